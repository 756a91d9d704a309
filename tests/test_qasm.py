"""OpenQASM 2.0 import (CPU): expressions, declarations, broadcasting, user
gates, errors, gate semantics against closed forms and brute force, and the
plans imported circuits get."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed, metrics, statevec as sv

qs = pytest.importorskip("paper_2609_19147_amd")
from paper_2609_19147_amd import qasm  # noqa: E402

HERE = os.path.join(os.path.dirname(__file__), "qasm")
HDR = 'OPENQASM 2.0;\ninclude "qelib1.inc";\n'


def as_oracle(gates):
    return [W.G(g.name, *g.wires, theta=g.theta, mat=g.mat) for g in gates]


def run(n, gates, psi0=None):
    psi0 = sv.basis(n, 0) if psi0 is None else psi0
    return sv.run(psi0, n, as_oracle(gates))


def one(src):
    n, g = qasm.loads(HDR + src)
    return n, g


@pytest.mark.parametrize("expr,val", [("pi/2", math.pi / 2), ("-pi/4", -math.pi / 4), ("2*pi/3", 2 * math.pi / 3),
                                      ("sin(pi/6)*2", 1.0), ("pi^2", math.pi ** 2), ("(1+2)*3", 9.0),
                                      ("1e-3", 1e-3), (".5", 0.5), ("-(-0.25)", 0.25), ("sqrt(4)+ln(exp(2))", 4.0),
                                      ("2^-1", 0.5), ("1-2-3", -4.0), ("8/2/2", 2.0)])
def test_expressions(expr, val):
    n, g = one(f"qreg q[1];\nrx({expr}) q[0];\n")
    assert g[0].name == "RX" and g[0].theta == pytest.approx(val, rel=1e-15, abs=1e-15)


def test_registers_broadcast_barrier_and_comments():
    n, g = one("qreg a[3];\nqreg b[3];\ncreg c[6];\n// comment\nh a;\nbarrier a,b;\ncx a, b;\ncz a[1], b;\n")
    assert n == 6
    assert [(x.name, x.wires) for x in g] == (
        [("H", (0,)), ("H", (1,)), ("H", (2,))] + [("CNOT", (k, 3 + k)) for k in range(3)]
        + [("CZ", (1, 3 + k)) for k in range(3)])


def test_files_load():
    n, g = qasm.load(os.path.join(HERE, "ghz_cat.qasm"), drop_measurements=True)
    assert n == 12 and sum(x.name == "CNOT" for x in g) == 10
    n, g = qasm.load(os.path.join(HERE, "user_gates.qasm"))
    assert n == 9 and len(g) > 30


@pytest.mark.parametrize("src,msg", [
    ("qreg q[2];\nfoo q[0];\n", "unknown gate"),
    ("qreg q[2];\ncx q[0];\n", "takes"),
    ("qreg q[2];\nrx q[0];\n", "takes"),
    ("qreg q[2];\ncx q[0], q[0];\n", "repeated"),
    ("qreg q[2];\nh q[2];\n", "out of range"),
    ("qreg q[2];\nh r[0];\n", "unknown register"),
    ("qreg q[2];\nqreg r[3];\ncx q, r;\n", "different sizes"),
    ("qreg q[2];\ncreg c[2];\nmeasure q -> c;\n", "not unitary"),
    ("qreg q[2];\nreset q[0];\n", "not unitary"),
    ("qreg q[2];\nopaque magic a;\nmagic q[0];\n", "opaque"),
    ("qreg q[2];\nrx(foo) q[0];\n", "unknown identifier"),
    ("qreg q[2];\nh q[0]\n", "missing ';'"),
])
def test_errors(src, msg):
    with pytest.raises(qasm.QasmError, match=msg):
        one(src)


def test_version_and_empty():
    with pytest.raises(qasm.QasmError):
        qasm.loads("OPENQASM 3.0;\nqreg q[1];\n")
    with pytest.raises(qasm.QasmError):
        qasm.loads(HDR)


def test_measurement_dropping():
    src = "qreg q[2];\ncreg c[2];\nh q[0];\ncx q[0],q[1];\nmeasure q -> c;\n"
    n, g = qasm.loads(HDR + src, drop_measurements=True)
    assert [x.name for x in g] == ["H", "CNOT"]
    with pytest.raises(qasm.QasmError, match="after a dropped measurement"):
        qasm.loads(HDR + src + "h q[1];\n", drop_measurements=True)


# ---------------------------------------------------------------- semantics
def mat_of(src, nq):
    """Full matrix of a small program by brute force over basis inputs."""
    n, g = one(f"qreg q[{nq}];\n" + src)
    cols = [run(n, g, sv.basis(n, j)) for j in range(1 << n)]
    return np.stack(cols, axis=1)


def test_single_qubit_definitions():
    th, ph, la = 0.7, -1.2, 0.4
    c, s = math.cos(th / 2), math.sin(th / 2)
    u3 = np.array([[c, -np.exp(1j * la) * s], [np.exp(1j * ph) * s, np.exp(1j * (ph + la)) * c]])
    assert np.allclose(mat_of(f"u3({th},{ph},{la}) q[0];\n", 1), u3, atol=1e-15)
    # u3(t, -pi/2, pi/2) = RX(t); u3(t, 0, 0) = RY(t); u2(f, l) = u3(pi/2, f, l); u1 = p = diag(1, e^il)
    assert np.allclose(mat_of(f"u3({th},-pi/2,pi/2) q[0];\n", 1), mat_of(f"rx({th}) q[0];\n", 1), atol=1e-15)
    assert np.allclose(mat_of(f"u3({th},0,0) q[0];\n", 1), mat_of(f"ry({th}) q[0];\n", 1), atol=1e-15)
    assert np.allclose(mat_of(f"u2({ph},{la}) q[0];\n", 1), mat_of(f"u3(pi/2,{ph},{la}) q[0];\n", 1), atol=1e-15)
    assert np.allclose(mat_of(f"u1({la}) q[0];\n", 1), np.diag([1, np.exp(1j * la)]), atol=1e-15)
    # rz differs from u1 by a global phase only
    rz, u1 = mat_of(f"rz({la}) q[0];\n", 1), mat_of(f"u1({la}) q[0];\n", 1)
    assert np.allclose(rz * np.exp(0.5j * la), u1, atol=1e-15)
    # sx^2 = x, sxdg sx = id
    assert np.allclose(mat_of("sx q[0];\nsx q[0];\n", 1), [[0, 1], [1, 0]], atol=1e-15)
    assert np.allclose(mat_of("sx q[0];\nsxdg q[0];\n", 1), np.eye(2), atol=1e-15)


def test_toffoli_and_fredkin_truth_tables():
    # qubit 0 is the most significant index bit
    T = mat_of("ccx q[0], q[1], q[2];\n", 3)
    F = mat_of("cswap q[0], q[1], q[2];\n", 3)
    for j in range(8):
        a, b, c = (j >> 2) & 1, (j >> 1) & 1, j & 1
        t = (a << 2) | (b << 1) | (c ^ (a & b))
        f = (a << 2) | ((c << 1) | b if a else (b << 1) | c)
        assert np.allclose(T[:, j], np.eye(8)[:, t], atol=1e-15)
        assert np.allclose(F[:, j], np.eye(8)[:, f], atol=1e-15)


def test_controlled_rotations():
    t = 0.9
    for name, U in (("crx", "rx"), ("cry", "ry"), ("crz", "rz")):
        M = mat_of(f"{name}({t}) q[0], q[1];\n", 2)
        u = mat_of(f"{U}({t}) q[0];\n", 1)
        assert np.allclose(M[:2, :2], np.eye(2), atol=1e-15) and np.allclose(M[2:, 2:], u, atol=1e-15)
        assert np.allclose(M[:2, 2:], 0) and np.allclose(M[2:, :2], 0)
    M = mat_of(f"cu1({t}) q[0], q[1];\n", 2)
    assert np.allclose(M, np.diag([1, 1, 1, np.exp(1j * t)]), atol=1e-15)


def qft_qasm(n):
    lines = [f"qreg q[{n}];"]
    for j in range(n):
        lines.append(f"h q[{j}];")
        for k in range(j + 1, n):
            lines.append(f"cu1(pi/{2 ** (k - j)}) q[{k}], q[{j}];")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("n", [3, 6, 9])
def test_qft_file_matches_closed_form(n):
    nq, g = one(qft_qasm(n))
    idx, c = W.sparse_state(n, 3, 4)
    psi0 = np.zeros(1 << n, complex)
    psi0[idx.astype(np.int64)] = c
    got = run(n, g, psi0)
    ref = closed.qft_sparse(n, idx, c, np.arange(1 << n, dtype=np.uint64))
    assert np.max(np.abs(got - ref)) < 1e-13


def test_ghz_file_state_and_plan():
    n, g = qasm.load(os.path.join(HERE, "ghz_cat.qasm"), drop_measurements=True)
    psi = run(n, g)
    # a: GHZ on qubits 0..6; b: cat state on qubits 7..11
    i0 = 0
    ia = sum(1 << (n - 1 - q) for q in range(7))
    ib = sum(1 << (n - 1 - q) for q in range(7, 12))
    ref = np.zeros(1 << n, complex)
    for x in (i0, ia, ib, ia | ib):
        ref[x] = 0.5
    assert np.max(np.abs(psi - ref)) < 1e-15
    # structured: each CNOT chain collapses into one permutation gather; the
    # default plan (dense windows allowed) needs no more layers than that
    kinds = [L["kind"] for L in qs.Plan(n, g, window_k=-1).describe()["layers"]]
    assert kinds.count("gf2") == 2 and "plain" not in kinds
    assert len(qs.Plan(n, g).describe()["layers"]) <= len(kinds)
    # one register alone: H pass + one gather
    src = "qreg q[10];\nh q[0];\n" + "".join(f"cx q[{k}],q[{k + 1}];\n" for k in range(9))
    n1, g1 = one(src)
    assert [L["kind"] for L in qs.Plan(n1, g1).describe()["layers"]] == ["tile", "gf2"]


def test_qft_file_fuses_like_the_native_stream():
    n = 16
    nq, g = one(qft_qasm(n))
    d = qs.Plan(n, g).describe()
    d0 = qs.Plan(n, W.qft_stream(n)).describe()
    assert [L["kind"] for L in d["layers"]] == [L["kind"] for L in d0["layers"]] == ["tile", "tile"]
    ops = [op["kind"] for L in d["layers"] for op in L["ops"]]
    assert ops == [op["kind"] for L in d0["layers"] for op in L["ops"]]


def test_user_gate_file_planned_exactly():
    from tests.plan_interp import run_plan
    n, g = qasm.load(os.path.join(HERE, "user_gates.qasm"))
    gates = as_oracle(g)
    psi0 = W.gaussian_state(n, 5)
    got = run_plan(qs.Plan(n, g).describe(), psi0, gates)
    assert np.max(np.abs(got - sv.run(psi0, n, gates))) < 1e-12
