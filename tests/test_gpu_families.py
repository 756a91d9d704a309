"""Weighted diagonal families on the GPU: long-range Ising Trotter steps (one
LUT group per bond distance) and the phase-estimation ladder with angles up
to 0.4 * 2^23 rad, against the oracle; the exact-phase QPE outcome at 21
qubits against its closed form."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import metrics, statevec as sv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


BAR = {"c64": 1e-10, "c128": 1e-24}


def run_both(qs, n, stream, dtype, psi0):
    st = qs.State(n, dtype, init=None)
    st.upload(psi0.astype(np.complex64 if dtype == "c64" else np.complex128))
    ref0 = st.download().astype(np.complex128)
    qs.apply(st, qs.Plan(n, stream))
    return st.download().astype(np.complex128), sv.run(ref0, n, stream)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_long_range_ising(qs, dtype):
    n = 12
    stream = W.long_range_ising_stream(n, 1.0, 1.5, 0.8, 0.05, 3)
    got, ref = run_both(qs, n, stream, dtype, W.gaussian_state(n, 4))
    assert metrics.infidelity(got, ref) <= BAR[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_qpe_ladder_large_angles(qs, dtype):
    t = 11
    stream = W.qpe_ladder_stream(t, 0.4, first_power=23 - (t - 1))
    got, ref = run_both(qs, t + 1, stream, dtype, sv.basis(t + 1, 0))
    assert metrics.infidelity(got, ref) <= BAR[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_qpe_exact_phase_21q(qs, dtype):
    t, j = 20, 704971
    st = qs.State(t + 1, dtype)
    qs.apply(st, qs.Plan(t + 1, W.qpe_ladder_stream(t, 2 * math.pi * j / 2 ** t)))
    amp = qs.amplitudes(st, [(j << 1) | 1])[0]
    assert abs(abs(amp) ** 2 - 1) < (1e-5 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_standalone_many_group_diagonal_layers(qs, dtype):
    """Diagonal-only streams become one standalone diagonal pass; with many
    groups it sums each amplitude's angle in FP64 (long-range ZZ couplings,
    13 distance groups; a controlled-power ladder with angles up to 0.4 2^23)."""
    n = 14
    lri = W.long_range_ising_stream(n, 1.0, 1.5, 0.0, 0.07, 1)[: n * (n - 1) // 2]
    ladder = [W.G("CPHASE", k, n - 1, theta=0.4 * 2.0 ** (10 + k)) for k in range(n - 1)]
    mixed = lri + ladder + [W.G("RZ", q, theta=0.3 + 0.1 * q) for q in range(n)]
    for stream in (lri, ladder, mixed):
        plan = qs.Plan(n, stream)
        assert [L["kind"] for L in plan.describe()["layers"]] == ["diag"]
        got, ref = run_both(qs, n, stream, dtype, W.gaussian_state(n, 6))
        assert metrics.infidelity(got, ref) <= BAR[dtype]
