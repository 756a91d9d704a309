"""XXZ / Heisenberg Trotter evolution and dense-window fusion on the GPU.

The open XXZ chain with a random field runs through the conjugated XX / YY
layers (one same-family run per Pauli pair); the two-leg ladder interleaves
XX, YY and ZZ per bond and runs as dense windows on the matrix cores; a QFT
written out as phase gates and CNOTs (no controlled-phase ladder left) and
random decomposed streams run as windows too.  All against the oracle at the
state bars (infidelity 1e-10 in complex64, 1e-24 in complex128); at 24 qubits
the window plan is checked against the structured plan of the same stream
and against the magnetisation the ladder conserves exactly.
"""
import numpy as np
import pytest

import workloads as W
from oracle import metrics, statevec as sv

pytestmark = pytest.mark.gpu

BAR = {"c64": 1e-10, "c128": 1e-24}


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


@pytest.fixture(autouse=True)
def _free_device_memory():
    yield
    import gc

    import torch
    gc.collect()
    torch.cuda.empty_cache()


def run_both(qs, n, stream, dtype, psi0, **opts):
    st = qs.State(n, dtype, init=None)
    st.upload(psi0.astype(np.complex64 if dtype == "c64" else np.complex128))
    ref0 = st.download().astype(np.complex128)
    plan = qs.Plan(n, stream, **opts)
    qs.apply(st, plan)
    return st, plan, st.download().astype(np.complex128), sv.run(ref0, n, stream), ref0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,delta", [(12, 1.0), (15, 0.5)])
def test_heisenberg_random_field_chain(qs, n, delta, dtype):
    stream = W.heisenberg_stream(n, 1.0, delta, 0.05, 3, W.random_fields(n, 1.0, n))
    st, plan, got, ref, _ = run_both(qs, n, stream, dtype, W.gaussian_state(n, 2))
    assert plan.describe()["windows"] == 0
    assert metrics.infidelity(got, ref) <= BAR[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("rungs,k", [(5, 0), (7, 4), (7, 6), (9, 5)])
def test_ladder_windows(qs, rungs, k, dtype):
    n = 2 * rungs
    stream = W.ladder_stream(rungs, 1.0, 0.5, 0.05, 2)
    st, plan, got, ref, psi0 = run_both(qs, n, stream, dtype, W.gaussian_state(n, rungs), window_k=k)
    d = plan.describe()
    assert d["windows"] > 0 and all(L["kind"] == "dense" for L in d["layers"])
    assert metrics.infidelity(got, ref) <= BAR[dtype]
    qs.apply(st, plan.inverse())
    assert metrics.infidelity(st.download().astype(np.complex128), psi0) <= BAR[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [10, 16])
def test_decomposed_qft(qs, n, dtype):
    stream = W.decomposed_qft_stream(n)
    st, plan, got, ref, _ = run_both(qs, n, stream, dtype, W.gaussian_state(n, 7))
    assert plan.describe()["windows"] > 0
    assert metrics.infidelity(got, ref) <= BAR[dtype]


@pytest.mark.parametrize("seed", range(4))
def test_random_decomposed_streams(qs, seed):
    n = 9 + seed
    stream = W.random_stream(n, 150, 70 + seed, kinds=("H", "RX", "RZ", "CNOT", "CZ", "SWAP", "RXX", "CU", "T"))
    for dtype in ("c64", "c128"):
        for k in (0, 4, 6):
            _, _, got, ref, _ = run_both(qs, n, stream, dtype, W.gaussian_state(n, seed), window_k=k)
            assert metrics.infidelity(got, ref) <= BAR[dtype], (dtype, k)


def test_ladder_24q_windows_match_structured_plan(qs):
    """24 qubits, one Trotter step from the Neel state: the dense-window plan
    and the structured plan (conjugated XX / YY layers in tile passes) agree,
    and both keep sum_q <Z_q> = 0 (each bond factor conserves it)."""
    rungs = 12
    n = 2 * rungs
    stream = W.ladder_stream(rungs, 1.0, 0.5, 0.05, 1)
    win = qs.Plan(n, stream)
    structured = qs.Plan(n, stream, window_k=-1)
    assert win.describe()["windows"] > 0 and structured.describe()["windows"] == 0
    a = qs.State(n, "c64")
    a.set_basis(W.neel_index(n))
    b = qs.State(n, "c64")
    b.set_basis(W.neel_index(n))
    qs.apply(a, win)
    qs.apply(b, structured)
    assert qs.infidelity(a, b) <= 1e-10
    for st in (a, b):
        assert abs(qs.expect(st, W.z_terms(n))) <= 1e-5
        assert abs(qs.norm2(st) - 1.0) <= 1e-5
