"""Imported OpenQASM 2.0 circuits on the GPU against the oracle (the same
gate list applied one gate at a time in complex128), at the state bars."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import metrics, statevec as sv

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(__file__), "qasm")
BAR = {"c64": 1e-10, "c128": 1e-24}


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


def check(qs, n, gates, dtype, **opts):
    psi0 = W.gaussian_state(n, 11).astype(np.complex64 if dtype == "c64" else np.complex128)
    st = qs.State(n, dtype, init=None)
    st.upload(psi0)
    qs.apply(st, qs.Plan(n, gates, **opts))
    ref = sv.run(psi0.astype(np.complex128), n, [W.G(g.name, *g.wires, theta=g.theta, mat=g.mat) for g in gates])
    assert metrics.infidelity(st.download().astype(np.complex128), ref) <= BAR[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("name", ["ghz_cat.qasm", "user_gates.qasm"])
@pytest.mark.parametrize("window_k", [0, -1])
def test_files(qs, name, dtype, window_k):
    from paper_2609_19147_amd import qasm
    n, g = qasm.load(os.path.join(HERE, name), drop_measurements=True)
    check(qs, n, g, dtype, window_k=window_k)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_qft_text_16q(qs, dtype):
    from paper_2609_19147_amd import qasm
    n = 16
    lines = ['OPENQASM 2.0;', 'include "qelib1.inc";', f"qreg q[{n}];"]
    for j in range(n):
        lines.append(f"h q[{j}];")
        lines += [f"cp(pi/{2 ** (k - j)}) q[{k}], q[{j}];" for k in range(j + 1, n)]
    nq, g = qasm.loads("\n".join(lines))
    check(qs, nq, g, dtype)
