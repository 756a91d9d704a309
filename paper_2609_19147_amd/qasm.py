"""OpenQASM 2.0 import (unitary subset).

The paper's import path reads OpenQASM 2.0 circuits, normalises gate names
into the detector vocabulary and skips barriers, so imported structured
circuits fuse as native ones do (Section "Benchmarks", QASM import, and
Appendix on the QASM sweep).  This reader covers the unitary part of the
language:

* ``OPENQASM 2.0;``, ``include "qelib1.inc";`` (the standard gates are
  built in), ``qreg`` (registers are numbered in declaration order), ``creg``;
* gate applications with parameter expressions (``pi``, ``+ - * / ^``, unary
  minus, ``sin cos tan exp ln sqrt``) and register broadcasting
  (``h q;``, ``cx a, b;`` over equal-size registers);
* user ``gate`` definitions, expanded on use; ``opaque`` declarations are
  rejected on use;
* ``barrier`` is skipped; ``measure``, ``reset`` and ``if`` are rejected
  (not unitary) unless ``drop_measurements`` is set, in which case trailing
  ``measure`` statements are dropped.

Gate names map onto the library's vocabulary: ``cx``/``CX`` -> CNOT,
``u1``/``p`` -> P, ``cu1``/``cp`` -> CPHASE, ``u2``/``u3``/``u``/``U`` -> U
(matrix), ``id`` -> I, controlled single-qubit gates -> CU (matrix of the
target block), ``ccx`` -> H, MCZ, H on the target, ``cswap`` -> CNOT, CCX,
CNOT.  ``rz`` is taken as exp(-i theta Z / 2) (qelib1's definition through
u1 differs by a global phase only).  Qubit q of the result is wire q of the
library (MSB-first: qubit 0 is the most significant index bit).
"""
from __future__ import annotations

import math
import re
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = ["QasmError", "QGate", "loads", "load"]


class QasmError(ValueError):
    pass


@dataclass(frozen=True)
class QGate:
    """One imported gate (the attributes the binding marshals)."""
    name: str
    wires: Tuple[int, ...]
    theta: float = 0.0
    param: int = -1
    scale: float = 1.0
    mat: Optional[Tuple[complex, ...]] = field(default=None, compare=False)

    def angle(self, params: Optional[Sequence[float]] = None) -> float:
        if self.param < 0:
            return float(self.theta)
        return float(self.theta) + float(self.scale) * float(params[self.param])


# ---------------------------------------------------------------- expressions
_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\.\d+(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)|([A-Za-z_]\w*)|(.))")
_FUNCS = {"sin": math.sin, "cos": math.cos, "tan": math.tan, "exp": math.exp, "ln": math.log, "sqrt": math.sqrt}


class _Expr:
    """Recursive-descent evaluator of OpenQASM 2.0 parameter expressions."""

    def __init__(self, text: str, env: Dict[str, float]):
        self.toks = []
        for num, name, op in _TOKEN.findall(text):
            if num:
                self.toks.append(("num", float(num)))
            elif name:
                self.toks.append(("name", name))
            elif op.strip():
                self.toks.append(("op", op))
        self.i = 0
        self.env = env

    def peek(self):
        return self.toks[self.i] if self.i < len(self.toks) else (None, None)

    def take(self, op=None):
        t = self.peek()
        if op is not None and t != ("op", op):
            raise QasmError(f"expected '{op}' in expression")
        self.i += 1
        return t

    def value(self) -> float:
        v = self.sum()
        if self.i != len(self.toks):
            raise QasmError("trailing tokens in expression")
        return v

    def sum(self) -> float:
        v = self.prod()
        while self.peek() in (("op", "+"), ("op", "-")):
            op = self.take()[1]
            r = self.prod()
            v = v + r if op == "+" else v - r
        return v

    def prod(self) -> float:
        v = self.unary()
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take()[1]
            r = self.unary()
            v = v * r if op == "*" else v / r
        return v

    def unary(self) -> float:
        if self.peek() == ("op", "-"):
            self.take()
            return -self.unary()
        if self.peek() == ("op", "+"):
            self.take()
            return self.unary()
        return self.power()

    def power(self) -> float:
        v = self.atom()
        if self.peek() == ("op", "^"):
            self.take()
            return v ** self.unary()
        return v

    def atom(self) -> float:
        kind, val = self.take()
        if kind == "num":
            return val
        if kind == "name":
            if val == "pi":
                return math.pi
            if val in _FUNCS:
                self.take("(")
                v = self.sum()
                self.take(")")
                return _FUNCS[val](v)
            if val in self.env:
                return self.env[val]
            raise QasmError(f"unknown identifier '{val}' in expression")
        if (kind, val) == ("op", "("):
            v = self.sum()
            self.take(")")
            return v
        raise QasmError("malformed expression")


def _split_top(text: str, sep: str = ",") -> List[str]:
    out, depth, cur = [], 0, []
    for ch in text:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == sep and depth == 0:
            out.append("".join(cur).strip())
            cur = []
        else:
            cur.append(ch)
    if "".join(cur).strip():
        out.append("".join(cur).strip())
    return out


# ---------------------------------------------------------------- matrices
def _u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]])


def _rx(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]])


def _ry(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -s], [s, c]])


def _rz(t):
    return np.diag([np.exp(-0.5j * t), np.exp(0.5j * t)])


_FIXED_1Q = {"h": np.array([[1, 1], [1, -1]]) / math.sqrt(2), "x": np.array([[0, 1], [1, 0]]),
             "y": np.array([[0, -1j], [1j, 0]]), "z": np.diag([1, -1]), "s": np.diag([1, 1j]),
             "sdg": np.diag([1, -1j]), "t": np.diag([1, np.exp(0.25j * math.pi)]),
             "tdg": np.diag([1, np.exp(-0.25j * math.pi)]),
             "sx": np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]]) / 2,
             "sxdg": np.array([[1 - 1j, 1 + 1j], [1 + 1j, 1 - 1j]]) / 2}


def _m(a: np.ndarray) -> Tuple[complex, ...]:
    return tuple(complex(v) for v in np.asarray(a, dtype=np.complex128).ravel())


# name -> (number of parameters, number of qubits)
_BUILTIN = {
    "id": (0, 1), "u0": (1, 1), "x": (0, 1), "y": (0, 1), "z": (0, 1), "h": (0, 1), "s": (0, 1),
    "sdg": (0, 1), "t": (0, 1), "tdg": (0, 1), "sx": (0, 1), "sxdg": (0, 1), "rx": (1, 1), "ry": (1, 1),
    "rz": (1, 1), "u1": (1, 1), "p": (1, 1), "u2": (2, 1), "u3": (3, 1), "u": (3, 1), "U": (3, 1),
    "cx": (0, 2), "CX": (0, 2), "cy": (0, 2), "cz": (0, 2), "ch": (0, 2), "csx": (0, 2), "swap": (0, 2),
    "crx": (1, 2), "cry": (1, 2), "crz": (1, 2), "cu1": (1, 2), "cp": (1, 2), "cu3": (3, 2), "cu": (4, 2),
    "rzz": (1, 2), "rxx": (1, 2), "ryy": (1, 2), "ccx": (0, 3), "cswap": (0, 3), "ccz": (0, 3),
}


def _builtin(name: str, p: Sequence[float], q: Sequence[int]) -> List[QGate]:
    if name == "id":
        return [QGate("I", (q[0],))]
    if name == "u0":
        return [QGate("I", (q[0],))]
    if name in ("x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx"):
        return [QGate(name.upper(), (q[0],))]
    if name == "sxdg":
        return [QGate("U", (q[0],), mat=_m(_FIXED_1Q["sxdg"]))]
    if name in ("rx", "ry", "rz"):
        return [QGate(name.upper(), (q[0],), theta=p[0])]
    if name in ("u1", "p"):
        return [QGate("P", (q[0],), theta=p[0])]
    if name == "u2":
        return [QGate("U", (q[0],), mat=_m(_u3(math.pi / 2, p[0], p[1])))]
    if name in ("u3", "u", "U"):
        return [QGate("U", (q[0],), mat=_m(_u3(p[0], p[1], p[2])))]
    if name in ("cx", "CX"):
        return [QGate("CNOT", (q[0], q[1]))]
    if name == "cz":
        return [QGate("CZ", (q[0], q[1]))]
    if name in ("cy", "ch", "csx"):
        return [QGate("CU", (q[0], q[1]), mat=_m(_FIXED_1Q[name[1:]]))]
    if name == "swap":
        return [QGate("SWAP", (q[0], q[1]))]
    if name in ("crx", "cry", "crz"):
        m = {"crx": _rx, "cry": _ry, "crz": _rz}[name](p[0])
        return [QGate("CU", (q[0], q[1]), mat=_m(m))]
    if name in ("cu1", "cp"):
        return [QGate("CPHASE", (q[0], q[1]), theta=p[0])]
    if name == "cu3":
        return [QGate("CU", (q[0], q[1]), mat=_m(_u3(p[0], p[1], p[2])))]
    if name == "cu":
        return [QGate("CU", (q[0], q[1]), mat=_m(np.exp(1j * p[3]) * _u3(p[0], p[1], p[2])))]
    if name in ("rzz", "rxx", "ryy"):
        return [QGate(name.upper(), (q[0], q[1]), theta=p[0])]
    if name == "ccz":
        return [QGate("MCZ", (q[0], q[1], q[2]))]
    if name == "ccx":
        return [QGate("H", (q[2],)), QGate("MCZ", (q[0], q[1], q[2])), QGate("H", (q[2],))]
    if name == "cswap":
        return ([QGate("CNOT", (q[2], q[1]))] + _builtin("ccx", (), (q[0], q[1], q[2]))
                + [QGate("CNOT", (q[2], q[1]))])
    raise QasmError(f"unknown gate '{name}'")


# ---------------------------------------------------------------- statements
@dataclass
class _GateDef:
    params: List[str]
    args: List[str]
    body: List[str]


_STMT_GATE = re.compile(r"^([A-Za-z_]\w*)\s*(?:\((.*)\))?\s+(.+)$", re.S)


def _strip_comments(text: str) -> str:
    return re.sub(r"//[^\n]*", "", text)


def _statements(text: str) -> List[str]:
    """Split into ';'-terminated statements, keeping gate bodies whole."""
    out, cur, depth = [], [], 0
    for ch in text:
        cur.append(ch)
        if ch == "{":
            depth += 1
        elif ch == "}":
            depth -= 1
            if depth == 0:
                out.append("".join(cur).strip())
                cur = []
        elif ch == ";" and depth == 0:
            out.append("".join(cur)[:-1].strip())
            cur = []
    if "".join(cur).strip():
        raise QasmError("missing ';' at the end of the program")
    return [s for s in out if s]


class _Reader:
    def __init__(self, drop_measurements: bool):
        self.regs: Dict[str, Tuple[int, int]] = {}
        self.nq = 0
        self.defs: Dict[str, _GateDef] = {}
        self.opaque = set()
        self.gates: List[QGate] = []
        self.drop_measurements = drop_measurements
        self.measured = False

    def operand(self, text: str) -> List[int]:
        m = re.fullmatch(r"\s*([A-Za-z_]\w*)\s*(?:\[\s*(\d+)\s*\])?\s*", text)
        if not m:
            raise QasmError(f"bad operand '{text}'")
        name, idx = m.group(1), m.group(2)
        if name not in self.regs:
            raise QasmError(f"unknown register '{name}'")
        off, size = self.regs[name]
        if idx is None:
            return list(range(off, off + size))
        if int(idx) >= size:
            raise QasmError(f"index {idx} out of range for '{name}'")
        return [off + int(idx)]

    def apply(self, name: str, params: List[float], qubits: List[int], depth: int = 0):
        if depth > 64:
            raise QasmError("gate definitions nest too deeply")
        if len(set(qubits)) != len(qubits):
            raise QasmError(f"repeated qubit in '{name}'")
        if name in self.defs:
            d = self.defs[name]
            if len(params) != len(d.params) or len(qubits) != len(d.args):
                raise QasmError(f"'{name}' takes {len(d.params)} parameters and {len(d.args)} qubits")
            env = dict(zip(d.params, params))
            amap = dict(zip(d.args, qubits))
            for st in d.body:
                nm, ps, ops = self.parse_app(st, env)
                sub = []
                for o in ops:
                    if o not in amap:
                        raise QasmError(f"unknown argument '{o}' in the body of '{name}'")
                    sub.append(amap[o])
                self.apply(nm, ps, sub, depth + 1)
            return
        if name in self.opaque:
            raise QasmError(f"opaque gate '{name}' has no definition")
        if name not in _BUILTIN:
            raise QasmError(f"unknown gate '{name}'")
        npar, nq = _BUILTIN[name]
        if len(params) != npar or len(qubits) != nq:
            raise QasmError(f"'{name}' takes {npar} parameters and {nq} qubits")
        self.gates.extend(_builtin(name, params, qubits))

    @staticmethod
    def parse_app(stmt: str, env: Dict[str, float]):
        m = _STMT_GATE.match(stmt.strip())
        if not m:
            raise QasmError(f"cannot parse '{stmt}'")
        name, ptext, otext = m.group(1), m.group(2), m.group(3)
        params = [_Expr(p, env).value() for p in _split_top(ptext)] if ptext and ptext.strip() else []
        ops = [o.strip() for o in otext.split(",")]
        return name, params, ops

    def statement(self, st: str):
        head = st.split(None, 1)[0] if st.split() else ""
        if st.startswith("OPENQASM"):
            if not re.fullmatch(r"OPENQASM\s+2(\.0)?", st):
                raise QasmError(f"unsupported version: '{st}'")
            return
        if head == "include":
            return  # the standard gates are built in
        if head in ("qreg", "creg"):
            m = re.fullmatch(r"(qreg|creg)\s+([A-Za-z_]\w*)\s*\[\s*(\d+)\s*\]", st)
            if not m:
                raise QasmError(f"bad declaration '{st}'")
            if m.group(1) == "qreg":
                if m.group(2) in self.regs:
                    raise QasmError(f"register '{m.group(2)}' declared twice")
                self.regs[m.group(2)] = (self.nq, int(m.group(3)))
                self.nq += int(m.group(3))
            return
        if head == "gate":
            m = re.fullmatch(r"gate\s+([A-Za-z_]\w*)\s*(?:\(([^)]*)\))?\s*([^{]*)\{(.*)\}", st, re.S)
            if not m:
                raise QasmError(f"bad gate definition '{st[:40]}'")
            params = [p.strip() for p in m.group(2).split(",")] if m.group(2) and m.group(2).strip() else []
            args = [a.strip() for a in m.group(3).split(",") if a.strip()]
            body = [b.strip() for b in m.group(4).split(";") if b.strip()]
            self.defs[m.group(1)] = _GateDef(params, args, [b for b in body if not b.startswith("barrier")])
            return
        if head == "opaque":
            m = re.match(r"opaque\s+([A-Za-z_]\w*)", st)
            self.opaque.add(m.group(1))
            return
        if head == "barrier":
            return
        if head == "measure":
            if self.drop_measurements:
                self.measured = True
                return
            raise QasmError("measure is not unitary (pass drop_measurements=True to drop trailing measurements)")
        if head in ("reset", "if"):
            raise QasmError(f"'{head}' is not unitary")
        if self.measured:
            raise QasmError("gate after a dropped measurement")
        name, params, ops = self.parse_app(st, {})
        regs = [self.operand(o) for o in ops]
        sizes = {len(r) for r in regs if len(r) > 1}
        if len(sizes) > 1:
            raise QasmError(f"registers of different sizes in '{st}'")
        width = sizes.pop() if sizes else 1
        for k in range(width):
            self.apply(name, params, [r[k] if len(r) > 1 else r[0] for r in regs])


def loads(text: str, drop_measurements: bool = False) -> Tuple[int, List[QGate]]:
    """Parse OpenQASM 2.0 source; returns (number of qubits, gates)."""
    R = _Reader(drop_measurements)
    for st in _statements(_strip_comments(text)):
        R.statement(" ".join(st.split()) if not st.startswith("gate") else st)
    if R.nq == 0:
        raise QasmError("no qubit register declared")
    return R.nq, R.gates


def load(path: str, drop_measurements: bool = False) -> Tuple[int, List[QGate]]:
    with open(path) as fh:
        return loads(fh.read(), drop_measurements)
