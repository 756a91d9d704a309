"""Dense k-qubit blocks (k = 4, 5, 6) on the matrix cores against the oracle.

Wire sets cover targets among the lowest state bits (the tile's column bits
then start above them), among the highest bits, interleaved, and random;
sizes span many tiles.  complex128 six-qubit blocks (matrix staged in LDS) are
checked the same way.  Bars as in the other parity tests.
"""
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


def run_device(qs, n, stream, dtype, seed=3):
    psi0 = W.gaussian_state(n, seed).astype(np.complex64 if dtype == "c64" else np.complex128)
    st = qs.State(n, dtype, init=None)
    st.upload(psi0)
    plan = qs.Plan(n, stream)
    qs.apply(st, plan)
    return st, plan, psi0.astype(np.complex128)


def check(got, ref, dtype, n):
    inf = metrics.infidelity(got, ref)
    assert inf <= (1e-10 if dtype == "c64" else 1e-24), inf
    amp = 1.0 / math.sqrt(1 << n)
    tol = (2e-5 if dtype == "c64" else 1e-12) * amp
    assert np.max(np.abs(got - ref)) <= tol, np.max(np.abs(got - ref)) / amp


def wire_sets(n, k):
    low = list(range(n - 1, n - 1 - k, -1))          # state bits 0..k-1
    high = list(range(k))                            # state bits n-k..n-1
    inter = list(range(0, 2 * k, 2))                 # every other bit from the top
    mixed = [n - 1, 0, n // 2, n - 3, 2, n // 2 + 1][:k]
    return [low, high, inter, mixed]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [4, 5, 6])
def test_structured_wire_sets(qs, k, dtype):
    n = 14
    rng = np.random.default_rng(100 + k)
    stream = [W.G("UNITARY", *w, mat=W.random_unitary(1 << k, rng)) for w in wire_sets(n, k)]
    st, plan, psi0 = run_device(qs, n, stream, dtype)
    assert [L["kind"] for L in plan.describe()["layers"]] == ["dense"] * 4
    check(st.download().astype(np.complex128), sv.run(psi0, n, stream), dtype, n)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k,n", [(4, 8), (4, 17), (5, 9), (5, 16), (6, 10), (6, 15)])
def test_random_blocks_with_other_layers(qs, k, n, dtype):
    stream = (W.dense_block_stream(n, 3, k, 7 * k + n) + W.qft_stream(n)
              + W.dense_block_stream(n, 2, k, 11 * k + n) + W.random_perm_block(n, 20, k))
    st, plan, psi0 = run_device(qs, n, stream, dtype)
    assert sum(L["kind"] == "dense" for L in plan.describe()["layers"]) == 5
    check(st.download().astype(np.complex128), sv.run(psi0, n, stream), dtype, n)
    # the inverse plan (conjugate-transposed blocks) returns the input
    qs.apply(st, plan.inverse())
    check(st.download().astype(np.complex128), psi0, dtype, n)


def test_dense_equals_plain_per_gate_path(qs):
    n, k = 16, 5
    stream = W.dense_block_stream(n, 6, k, 77)
    st, plan, psi0 = run_device(qs, n, stream, "c64")
    ref = qs.State(n, "c64", init=None)
    ref.upload(psi0.astype(np.complex64))
    qs.apply_gates(ref, stream)
    assert qs.infidelity(st, ref) <= 1e-10


@pytest.mark.parametrize("dtype,k", [("c64", 6), ("c64", 5), ("c128", 6)])
def test_many_tile_blocks_at_24_qubits_against_oracle(qs, dtype, k):
    """24 qubits (2^18 tiles over the persistent grid, each workgroup walking
    a hundred tiles, as at the benchmark's 30 qubits): three seeded k-qubit
    blocks against the oracle, element by element, then the inverse plan
    back to the input and the norm."""
    n = 24
    stream = W.dense_block_stream(n, 3, k, 500 + k)
    st, plan, psi0 = run_device(qs, n, stream, dtype, seed=9)
    assert [L["kind"] for L in plan.describe()["layers"]] == ["dense"] * 3
    check(st.download().astype(np.complex128), sv.run(psi0, n, stream), dtype, n)
    qs.apply(st, plan.inverse())
    check(st.download().astype(np.complex128), psi0, dtype, n)
    assert abs(qs.norm2(st) - metrics.norm2(psi0)) <= (1e-6 if dtype == "c64" else 1e-13)
