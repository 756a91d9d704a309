"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* inputs: gate streams (lists of :class:`Gate`),
Pauli observables (lists of ``(coeff, x_mask, z_mask)``), graphs and seeded
random states.  It contains none of the simulation arithmetic: it never
applies a gate, never forms a matrix product and never evaluates an
expectation.  Both the CPU oracle (``oracle/``) and the HIP path
(``paper_2609_19147_amd``) consume exactly what is produced here.

Conventions (Section "State Management" and the gate-operation description
of the paper): qubit ``q`` is bit ``n-1-q`` of the basis index (MSB-first).
Pauli masks use *qubit* numbering: bit ``q`` of ``x_mask``/``z_mask`` refers
to qubit ``q``; a qubit with both bits set carries a Y.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate names understood by both sides.  Matrices are defined by the oracle
# (the plain definition) and independently by the library.
ONE_QUBIT = ("I", "H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX",
             "RX", "RY", "RZ", "P", "U")
TWO_QUBIT = ("CNOT", "CZ", "CPHASE", "SWAP", "RZZ", "RXX", "RYY", "CU")
MULTI = ("MCZ", "MCP", "UNITARY")
PARAMETRIC = ("RX", "RY", "RZ", "P", "CPHASE", "RZZ", "RXX", "RYY", "MCP")


@dataclass(frozen=True)
class Gate:
    """One gate of a stream.

    ``wires`` lists qubits (for controlled gates: control(s) first, target
    last).  ``theta`` is the fixed angle.  When ``param >= 0`` the angle is
    ``theta + scale * params[param]`` (parameters are bound at run time).
    ``mat`` is a row-major complex matrix for ``U`` (2x2), ``CU`` (the
    2x2 target block) and ``UNITARY`` (2^k x 2^k, first wire = most
    significant row bit).
    """
    name: str
    wires: Tuple[int, ...]
    theta: float = 0.0
    param: int = -1
    scale: float = 1.0
    mat: Optional[Tuple[complex, ...]] = field(default=None, compare=False)

    def angle(self, params: Optional[Sequence[float]] = None) -> float:
        if self.param < 0:
            return float(self.theta)
        if params is None:
            raise ValueError(f"gate {self.name} needs parameter {self.param}")
        return float(self.theta) + float(self.scale) * float(params[self.param])


def G(name: str, *wires: int, theta: float = 0.0, param: int = -1,
      scale: float = 1.0, mat=None) -> Gate:
    m = None if mat is None else tuple(complex(v) for v in np.asarray(mat).ravel())
    return Gate(name, tuple(int(w) for w in wires), float(theta), int(param),
                float(scale), m)


# --------------------------------------------------------------------------
# Seeded states
# --------------------------------------------------------------------------

def gaussian_state(n: int, seed: int) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes, normalised in FP64 (complex128).

    ``numpy.random.default_rng(seed)`` (PCG64); real parts are drawn first,
    then imaginary parts.  Callers that run in complex64 cast this array and
    hand the *rounded* values (upcast) to the oracle.
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(1 << n)
    im = rng.standard_normal(1 << n)
    psi = re + 1j * im
    psi /= math.sqrt(float(np.vdot(psi, psi).real))
    return psi


def sparse_state(n: int, seed: int, k: int = 8) -> Tuple[np.ndarray, np.ndarray]:
    """``k`` distinct random basis indices with random complex weights.

    Returns ``(indices, coeffs)`` (uint64, complex128), coefficients
    normalised.  Used at sizes where a dense host state is too large: every
    output amplitude of a linear map is then a ``k``-term sum.
    """
    rng = np.random.default_rng(seed)
    idx = np.unique(rng.integers(0, 1 << n, size=4 * k, dtype=np.uint64))[:k]
    rng.shuffle(idx)
    c = rng.standard_normal(len(idx)) + 1j * rng.standard_normal(len(idx))
    c /= math.sqrt(float(np.vdot(c, c).real))
    return idx.astype(np.uint64), c


def index_tag_state(n: int) -> np.ndarray:
    """State whose amplitude at index i encodes i exactly in complex64.

    Re = i mod 2^24, Im = floor(i / 2^24); both are integers below 2^24 and
    therefore exact in float32.  Not normalised: it is a probe for
    permutations, which move amplitudes without arithmetic.
    """
    i = np.arange(1 << n, dtype=np.int64)
    return ((i & ((1 << 24) - 1)).astype(np.float64)
            + 1j * (i >> 24).astype(np.float64))


# --------------------------------------------------------------------------
# Gate streams
# --------------------------------------------------------------------------

def qft_stream(n: int) -> List[Gate]:
    """Textbook QFT: for j: H(j), then CPHASE(pi/2^(k-j)) on (k, j), k>j.

    No final swaps, so the output is bit-reversed; n + n(n-1)/2 gates
    (Section "Quantum Fourier Transform" and the benchmark depth formulas).
    """
    out: List[Gate] = []
    for j in range(n):
        out.append(G("H", j))
        for k in range(j + 1, n):
            out.append(G("CPHASE", k, j, theta=math.pi / (1 << (k - j))))
    return out


def qft_register_stream(qubits: Sequence[int], degree: Optional[int] = None) -> List[Gate]:
    """QFT stream on the listed qubits (most significant first), no swaps.

    Same gate order as :func:`qft_stream`, with register position ``j``
    standing for ``qubits[j]``.  ``degree`` keeps only the controlled phases
    whose register distance ``k - j`` is at most ``degree`` (the approximate
    QFT); ``None`` keeps them all.
    """
    out: List[Gate] = []
    m = len(qubits)
    for j in range(m):
        out.append(G("H", qubits[j]))
        for k in range(j + 1, m):
            if degree is not None and k - j > degree:
                break
            out.append(G("CPHASE", qubits[k], qubits[j], theta=math.pi / (1 << (k - j))))
    return out


def wht_stream(n: int) -> List[Gate]:
    return [G("H", q) for q in range(n)]


def random_perm_block(n: int, n_gates: int, seed: int) -> List[Gate]:
    """Random X / CNOT / SWAP block: kind uniform, wires uniform distinct."""
    rng = np.random.default_rng(seed)
    out: List[Gate] = []
    for _ in range(n_gates):
        kind = int(rng.integers(0, 3))
        w = rng.choice(n, size=2, replace=False)
        if kind == 0:
            out.append(G("X", int(w[0])))
        elif kind == 1:
            out.append(G("CNOT", int(w[0]), int(w[1])))
        else:
            out.append(G("SWAP", int(w[0]), int(w[1])))
    return out


def ghz_stream(n: int) -> List[Gate]:
    return [G("H", 0)] + [G("CNOT", q, q + 1) for q in range(n - 1)]


def tfim_first_order_stream(n: int, J: float, h: float, t: float, r: int) -> List[Gate]:
    """First-order Lie-Trotter TFIM (open chain), ZZ layer before X layer.

    H = -J sum Z_i Z_{i+1} + h sum X_i; exp(i J Z Z dt) = RZZ(-2 J dt) and
    exp(-i h X dt) = RX(2 h dt), dt = t / r; start |0...0>.
    """
    dt = t / r
    out: List[Gate] = []
    for _ in range(r):
        out += [G("RZZ", q, q + 1, theta=-2.0 * J * dt) for q in range(n - 1)]
        out += [G("RX", q, theta=2.0 * h * dt) for q in range(n)]
    return out


def tfim_strang_stream(n: int, J: float, h: float, dt: float, steps: int,
                       h_layer: bool = True) -> List[Gate]:
    """Second-order (Strang) TFIM steps: RX(h dt), RZZ(-2 J dt), RX(h dt).

    Optionally preceded by an H layer on every qubit.
    """
    out: List[Gate] = wht_stream(n) if h_layer else []
    for _ in range(steps):
        out += [G("RX", q, theta=h * dt) for q in range(n)]
        out += [G("RZZ", q, q + 1, theta=-2.0 * J * dt) for q in range(n - 1)]
        out += [G("RX", q, theta=h * dt) for q in range(n)]
    return out


def hea_stream(n: int, layers: int) -> List[Gate]:
    """Hardware-efficient ansatz: per layer RY then RZ on every qubit, then
    CNOT(q, q+1) for q = 0..n-2.  Parameter index = (layer*n + q)*2 + {0: RY, 1: RZ}.
    """
    out: List[Gate] = []
    for l in range(layers):
        for q in range(n):
            out.append(G("RY", q, param=(l * n + q) * 2))
            out.append(G("RZ", q, param=(l * n + q) * 2 + 1))
        out += [G("CNOT", q, q + 1) for q in range(n - 1)]
    return out


def hea_params(n: int, layers: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-math.pi, math.pi, size=2 * n * layers)


def random_regular3_graph(n: int, rng: np.random.Generator) -> List[Tuple[int, int]]:
    """Random 3-regular simple graph: configuration model with rejection."""
    if (3 * n) % 2:
        raise ValueError("a 3-regular graph needs an even vertex count")
    while True:
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted(seen)


@dataclass
class QaoaInstance:
    n: int
    edges: List[Tuple[int, int]]
    gammas: np.ndarray
    betas: np.ndarray


def qaoa_instances(count: int, seed: int, depth: int = 4,
                   n_choices: Sequence[int] = (16, 18, 20, 22, 24)) -> List[QaoaInstance]:
    """MaxCut QAOA instances: n uniform over ``n_choices`` (even, so that a
    3-regular graph exists), random 3-regular graph, gamma, beta ~ U[0, pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(n_choices)))
        edges = random_regular3_graph(n, rng)
        gam = rng.uniform(0.0, math.pi, size=depth)
        bet = rng.uniform(0.0, math.pi, size=depth)
        out.append(QaoaInstance(n, edges, gam, bet))
    return out


def qaoa_stream(inst: QaoaInstance, param_offset: int = -1, h_layer: bool = True) -> List[Gate]:
    """|+>^n (an H layer on |0...0>, omitted with ``h_layer=False`` for runs
    that start from |+>^n directly), then per layer exp(-i gamma C) (as
    RZZ(-gamma) per edge, equal to the cost unitary up to a global phase) and
    exp(-i beta sum X) = RX(2 beta).

    With ``param_offset >= 0`` the angles are parameters: gamma_l at index
    offset + 2l (RZZ scale -1), beta_l at offset + 2l + 1 (RX scale 2).
    """
    out = wht_stream(inst.n) if h_layer else []
    for l in range(len(inst.gammas)):
        if param_offset >= 0:
            out += [G("RZZ", u, v, param=param_offset + 2 * l, scale=-1.0) for u, v in inst.edges]
            out += [G("RX", q, param=param_offset + 2 * l + 1, scale=2.0) for q in range(inst.n)]
        else:
            out += [G("RZZ", u, v, theta=-float(inst.gammas[l])) for u, v in inst.edges]
            out += [G("RX", q, theta=2.0 * float(inst.betas[l])) for q in range(inst.n)]
    return out


def grover_stream(n: int, marked: int, iterations: int) -> List[Gate]:
    """Grover search: H layer, then per iteration an oracle (X-conjugated
    multi-controlled Z marking ``marked``, given MSB-first) and the diffusion
    H X MCZ X H."""
    allq = tuple(range(n))
    zeros = [q for q in range(n) if not (marked >> (n - 1 - q)) & 1]
    out = wht_stream(n)
    for _ in range(iterations):
        out += [G("X", q) for q in zeros]
        out.append(G("MCZ", *allq))
        out += [G("X", q) for q in zeros]
        out += wht_stream(n)
        out += [G("X", q) for q in range(n)]
        out.append(G("MCZ", *allq))
        out += [G("X", q) for q in range(n)]
        out += wht_stream(n)
    return out


# --------------------------------------------------------------------------
# Observables: lists of (coeff, x_mask, z_mask), bit q = qubit q
# --------------------------------------------------------------------------

PauliTerm = Tuple[float, int, int]


def pauli(coeff: float, ops: dict) -> PauliTerm:
    """``ops`` maps qubit -> 'X' | 'Y' | 'Z'."""
    xm = zm = 0
    for q, p in ops.items():
        if p in ("X", "Y"):
            xm |= 1 << q
        if p in ("Z", "Y"):
            zm |= 1 << q
    return (float(coeff), xm, zm)


def xxz_terms(n: int, jz: float = 0.5, J: float = 1.0) -> List[PauliTerm]:
    """Open-chain XXZ: J sum_i (X_i X_{i+1} + Y_i Y_{i+1} + jz Z_i Z_{i+1})."""
    out: List[PauliTerm] = []
    for i in range(n - 1):
        out.append(pauli(J, {i: "X", i + 1: "X"}))
        out.append(pauli(J, {i: "Y", i + 1: "Y"}))
        out.append(pauli(J * jz, {i: "Z", i + 1: "Z"}))
    return out


def z_terms(n: int) -> List[PauliTerm]:
    return [pauli(1.0, {q: "Z"}) for q in range(n)]


def x_terms(n: int) -> List[PauliTerm]:
    return [pauli(1.0, {q: "X"}) for q in range(n)]


def zz_chain_terms(n: int) -> List[PauliTerm]:
    return [pauli(1.0, {q: "Z", q + 1: "Z"}) for q in range(n - 1)]


def maxcut_terms(edges: Sequence[Tuple[int, int]]) -> List[PauliTerm]:
    """C = sum_E (1 - Z_u Z_v) / 2 as Pauli terms (identity term has masks 0)."""
    out: List[PauliTerm] = [(0.5 * len(edges), 0, 0)]
    out += [pauli(-0.5, {u: "Z", v: "Z"}) for u, v in edges]
    return out


def random_stream(n: int, n_gates: int, seed: int, kinds: Sequence[str] = None) -> List[Gate]:
    """Random mixed stream over the whole vocabulary (for parity tests)."""
    rng = np.random.default_rng(seed)
    kinds = list(kinds or ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY",
                           "RZ", "P", "U", "CNOT", "CZ", "CPHASE", "SWAP", "RZZ", "RXX",
                           "RYY", "CU"))
    out: List[Gate] = []
    for _ in range(n_gates):
        k = kinds[int(rng.integers(0, len(kinds)))]
        th = float(rng.uniform(-math.pi, math.pi))
        if k in ONE_QUBIT:
            q = int(rng.integers(0, n))
            if k == "U":
                out.append(G("U", q, mat=random_unitary(2, rng)))
            else:
                out.append(G(k, q, theta=th))
        else:
            w = rng.choice(n, size=2, replace=False)
            if k == "CU":
                out.append(G("CU", int(w[0]), int(w[1]), mat=random_unitary(2, rng)))
            else:
                out.append(G(k, int(w[0]), int(w[1]), theta=th))
    return out


def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-ish unitary: QR of a complex Gaussian matrix, phases fixed.

    (Input generation only: the result is a list of numbers handed to both
    sides as a gate matrix.)"""
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))


def long_range_ising_stream(n: int, j0: float, alpha: float, h: float, dt: float, steps: int) -> List[Gate]:
    """Long-range transverse-field Ising Trotter evolution from |0...0>:
    H = -sum_{i<j} J(|i-j|) Z_i Z_j + h sum_i X_i with J(r) = j0 / r^alpha (all
    n(n-1)/2 bonds, n-1 distance classes).  Per first-order step: the ZZ layer
    as RZZ(-2 J(r) dt) on every bond (bonds ordered by distance), then
    RX(2 h dt) on every qubit."""
    out: List[Gate] = []
    for _ in range(steps):
        for r in range(1, n):
            th = -2.0 * j0 / r ** alpha * dt
            out += [G("RZZ", i, i + r, theta=th) for i in range(n - r)]
        out += [G("RX", q, theta=2.0 * h * dt) for q in range(n)]
    return out


def qpe_ladder_stream(t: int, theta: float, first_power: int = 0) -> List[Gate]:
    """Phase estimation of P(theta) on one target qubit (wire t, prepared in
    |1>, its e^{i theta} eigenstate) with t counting qubits: H on the counting
    wires, controlled-P(theta 2^(first_power + k)) from counting wire k to the
    target, then the inverse QFT (the QFT stream reversed, conjugated) on the
    counting wires.  For theta 2^first_power = 2 pi j / 2^t the counting
    register ends in |j> exactly.  The ladder's angles reach
    theta 2^(first_power + t - 1)."""
    out: List[Gate] = [G("X", t)] + [G("H", q) for q in range(t)]
    for k in range(t):
        out.append(G("CPHASE", k, t, theta=theta * 2.0 ** (first_power + k)))
    inv = []
    for g in reversed(qft_stream(t)):
        inv.append(G("CPHASE", *g.wires, theta=-g.theta) if g.name == "CPHASE" else g)
    return out + inv


def random_fields(n: int, width: float, seed: int) -> np.ndarray:
    """Random longitudinal fields h_q ~ U[-width, width] (seeded)."""
    return np.random.default_rng(seed).uniform(-width, width, size=n)


def heisenberg_stream(n: int, J: float, delta: float, dt: float, steps: int,
                      fields: Optional[Sequence[float]] = None) -> List[Gate]:
    """First-order Trotter evolution under the open-chain XXZ Hamiltonian
    H = J sum_i (X_i X_{i+1} + Y_i Y_{i+1} + delta Z_i Z_{i+1}) + sum_q h_q Z_q.
    Per step: RXX(2 J dt) on every bond, then RYY(2 J dt) on every bond, then
    RZZ(2 J delta dt) on every bond, then RZ(2 h_q dt) per qubit (one same-family
    run per Pauli pair; delta = 1 is the Heisenberg chain)."""
    out: List[Gate] = []
    for _ in range(steps):
        for name, th in (("RXX", 2.0 * J * dt), ("RYY", 2.0 * J * dt), ("RZZ", 2.0 * J * delta * dt)):
            out += [G(name, i, i + 1, theta=th) for i in range(n - 1)]
        if fields is not None:
            out += [G("RZ", q, theta=2.0 * float(fields[q]) * dt) for q in range(n)]
    return out


def ladder_bonds(rungs: int) -> List[Tuple[int, int]]:
    """Bonds of a two-leg ladder with site (rung r, leg l) on qubit 2 r + l, in
    rung order: the rung (2r, 2r+1), then the leg bonds to rung r + 1."""
    out: List[Tuple[int, int]] = []
    for r in range(rungs):
        out.append((2 * r, 2 * r + 1))
        if r + 1 < rungs:
            out += [(2 * r, 2 * r + 2), (2 * r + 1, 2 * r + 3)]
    return out


def ladder_stream(rungs: int, J: float, delta: float, dt: float, steps: int) -> List[Gate]:
    """First-order Trotter evolution of the two-leg XXZ ladder
    H = J sum_bonds (XX + YY + delta ZZ): per step and per bond, in bond order,
    RXX(2 J dt), RYY(2 J dt), RZZ(2 J delta dt).  The three Pauli pairs of one
    bond commute, so each bond's triple is exactly exp(-i dt h_bond); the
    families interleave, so no same-family run forms."""
    out: List[Gate] = []
    for _ in range(steps):
        for a, b in ladder_bonds(rungs):
            out += [G("RXX", a, b, theta=2.0 * J * dt), G("RYY", a, b, theta=2.0 * J * dt),
                    G("RZZ", a, b, theta=2.0 * J * delta * dt)]
    return out


def neel_index(n: int) -> int:
    """Basis index of |0101...> (qubit q in state q mod 2)."""
    return sum(1 << (n - 1 - q) for q in range(1, n, 2))


def decomposed_qft_stream(n: int) -> List[Gate]:
    """The QFT stream with every controlled phase written out as phase gates
    and CNOTs: CP(t) on (c, g) = P(t/2) c, CNOT(c, g), P(-t/2) g, CNOT(c, g),
    P(t/2) g (the form a transpiled file carries; no controlled-phase ladder
    remains for a stage detector)."""
    out: List[Gate] = []
    for g in qft_stream(n):
        if g.name != "CPHASE":
            out.append(g)
            continue
        c, t = g.wires
        th = g.theta
        out += [G("P", c, theta=th / 2), G("CNOT", c, t), G("P", t, theta=-th / 2), G("CNOT", c, t),
                G("P", t, theta=th / 2)]
    return out


def dense_block_stream(n: int, count: int, k: int, seed: int) -> List[Gate]:
    """``count`` UNITARY gates on k distinct random wires each, with Haar-ish
    2^k x 2^k matrices (the dense-block microbenchmark's input)."""
    rng = np.random.default_rng(seed)
    out: List[Gate] = []
    for _ in range(count):
        w = rng.choice(n, size=k, replace=False)
        out.append(G("UNITARY", *[int(x) for x in w], mat=random_unitary(1 << k, rng)))
    return out


def gaussian_state_torch(n: int, seed: int, dtype: str = "c64", out=None):
    """Seeded i.i.d. complex Gaussian state generated on the GPU with torch's
    Philox generator, normalised in FP64 (for sizes where a host state would be
    impractical, e.g. 30 qubits).  Writes into ``out`` when given."""
    import torch
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    psi = out if out is not None else torch.empty(1 << n, dtype=tdt, device="cuda")
    chunk = 1 << 26
    for s in range(0, 1 << n, chunk):
        psi[s:s + chunk] = torch.randn(min(chunk, (1 << n) - s), dtype=tdt, device="cuda", generator=g)
    nrm = torch.linalg.vector_norm(psi.view(torch.float32 if dtype == "c64" else torch.float64), dtype=torch.float64)
    psi /= nrm.to(psi.real.dtype)
    return psi
