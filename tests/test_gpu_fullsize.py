"""Full-size parity: the state-vector benchmark's circuit and launch
configuration at 30 qubits, the 25-qubit TFIM evolution, and a 30-qubit GF(2)
permutation, checked on sampled outputs that the oracle computes one by one
(closed forms, a stored oracle run) and on properties that hold at any size.

Bars: relative L2 error over the sampled amplitudes <= 1e-5 in complex64 and
<= 1e-12 in complex128 (the square roots of the infidelity bars 1e-10 and
1e-24); permutations bit-exact.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REL = {"c64": 1e-5, "c128": 1e-12}
N30 = 30


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


def rel_err(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def sparse_on_device(qs, n, dtype, seed, k=8):
    """A k-sparse state written straight into device memory; returns the
    coefficients as the device holds them (rounded to the dtype)."""
    import torch
    idx, c = W.sparse_state(n, seed, k)
    nd = np.complex64 if dtype == "c64" else np.complex128
    c = c.astype(nd)
    st = qs.State(n, dtype, init=None)
    t = st.tensor()
    t.zero_()
    t[torch.as_tensor(idx.astype(np.int64), device="cuda")] = torch.as_tensor(c, device="cuda")
    return st, idx, c.astype(np.complex128)


def sample_indices(n, seed, count=8192):
    rng = np.random.default_rng(seed)
    ys = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return np.unique(np.concatenate([ys, np.array([0, (1 << n) - 1], np.uint64)]))


@pytest.mark.parametrize("dtype,tile_bits", [("c64", 0), ("c128", 0), ("c64", 14), ("c128", 12), ("c64", 12)])
def test_benchmark_circuit_30q_sampled_outputs(qs, dtype, tile_bits):
    """The benchmark's plan (same circuit, same planner options) on a sparse
    input: out[y] = (Walsh . QFT psi0)[src(y)] with src from the X/CNOT/SWAP block.
    Tiles that fill the LDS (2^13 complex128, 2^14 complex64 amplitudes) run
    the pipelined kernel, one workgroup per CU walking 512 cosets."""
    from bench import BLOCK_SEED, circuit
    stream = circuit(N30)
    plan = qs.Plan(N30, stream, max_tile_bits=tile_bits)
    kinds = [L["kind"] for L in plan.describe()["layers"]]
    assert kinds[-1] == "gf2" and set(kinds[:-1]) == {"tile"}
    assert len(kinds) == (5 if tile_bits == 12 else 4)
    st, idx, c = sparse_on_device(qs, N30, dtype, seed=5)
    qs.apply(st, plan)
    ys = sample_indices(N30, 11)
    got = qs.amplitudes(st, ys).astype(np.complex128)
    perm = W.random_perm_block(N30, 200, BLOCK_SEED)
    assert stream[-200:] == perm
    ref = closed.qft_wht_sparse(N30, idx, c, closed.perm_source(N30, perm, ys))
    assert rel_err(got, ref) <= REL[dtype], rel_err(got, ref)
    # the whole state keeps its norm
    assert abs(qs.norm2(st) - float(np.vdot(c, c).real)) <= (1e-5 if dtype == "c64" else 1e-12)


def test_benchmark_input_round_trip_30q(qs):
    """The benchmark's exact input (seeded Gaussian, 30 qubits, complex64):
    the plan followed by its inverse plan returns it."""
    from bench import STATE_SEED, circuit
    plan = qs.Plan(N30, circuit(N30))
    st = qs.State(N30, "c64", init=None)
    W.gaussian_state_torch(N30, STATE_SEED, "c64", out=st.tensor())
    ref = qs.State(N30, "c64", init=None, lazy_scratch=True)
    ref.copy_from(st)
    n0 = qs.norm2(st)
    qs.apply(st, plan)
    assert abs(qs.norm2(st) - n0) <= 1e-5
    qs.apply(st, plan.inverse())
    assert qs.infidelity(st, ref) <= 1e-10


def test_gf2_block_30q_index_tags_bit_exact(qs):
    """The benchmark's 200-gate X/CNOT/SWAP block as one GF(2) gather at 30
    qubits on a state whose amplitude at i encodes i exactly."""
    import torch
    from bench import BLOCK_SEED
    perm = W.random_perm_block(N30, 200, BLOCK_SEED)
    plan = qs.Plan(N30, perm)
    assert [L["kind"] for L in plan.describe()["layers"]] == ["gf2"]
    st = qs.State(N30, "c64", init=None)
    t = st.tensor()
    chunk = 1 << 26
    for s in range(0, 1 << N30, chunk):
        i = torch.arange(s, s + chunk, dtype=torch.int64, device="cuda")
        t[s:s + chunk] = torch.complex((i & ((1 << 24) - 1)).to(torch.float32), (i >> 24).to(torch.float32))
    qs.apply(st, plan)
    ys = sample_indices(N30, 17, 65536)
    got = qs.amplitudes(st, ys)
    src = closed.perm_source(N30, perm, ys)
    want = ((src & np.uint64((1 << 24) - 1)).astype(np.float32)
            + 1j * (src >> np.uint64(24)).astype(np.float32)).astype(np.complex64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_tfim25_strang_against_stored_oracle_run(qs, dtype):
    """25-qubit open-chain TFIM (J = 1, h = 0.8, dt = 0.05, 40 Strang steps from
    the H layer on |0...0>) against the oracle's stored run: sampled amplitudes,
    <X_i>, <Z_i Z_i+1>, and <Z_i> = 0 (the global spin flip commutes with H and
    fixes the initial state)."""
    with open(os.path.join(HERE, "golden", "tfim25_strang.json")) as fh:
        gold = json.load(fh)
    w = gold["workload"]
    stream = W.tfim_strang_stream(w["n"], w["J"], w["h"], w["dt"], w["steps"])
    assert len(stream) == w["gates"]
    plan = qs.Plan(w["n"], stream)
    st = qs.State(w["n"], dtype)
    qs.apply(st, plan)
    got = qs.amplitudes(st, np.array(gold["sample_idx"], np.uint64)).astype(np.complex128)
    ref = np.array(gold["sample_re"]) + 1j * np.array(gold["sample_im"])
    assert rel_err(got, ref) <= REL[dtype], rel_err(got, ref)
    obs_tol = 2e-5 if dtype == "c64" else 1e-11
    _, x = qs.expect(st, W.x_terms(w["n"]), per_term=True)
    _, zz = qs.expect(st, W.zz_chain_terms(w["n"]), per_term=True)
    _, z = qs.expect(st, W.z_terms(w["n"]), per_term=True)
    assert np.max(np.abs(x - np.array(gold["x"]))) <= obs_tol
    assert np.max(np.abs(zz - np.array(gold["zz"]))) <= obs_tol
    assert np.max(np.abs(z)) <= obs_tol
    assert abs(qs.norm2(st) - 1.0) <= (1e-5 if dtype == "c64" else 1e-12)


def test_max_qubits_32_benchmark_shape(qs):
    """The largest state the library takes (32 qubits, 32 GiB complex64 plus an
    equal gather buffer): QFT -> Walsh -> 60-gate X/CNOT/SWAP block on a sparse
    input, sampled outputs against the closed form, the norm fused into the
    gather, and the block alone on index tags bit for bit."""
    import torch
    n = 32
    perm = W.random_perm_block(n, 60, 33)
    stream = W.qft_stream(n) + W.wht_stream(n) + perm
    plan = qs.Plan(n, stream)
    assert [L["kind"] for L in plan.describe()["layers"]][-1] == "gf2"
    st, idx, c = sparse_on_device(qs, n, "c64", seed=9)
    nrm = qs.apply_norm2(st, plan)
    assert abs(nrm - float(np.vdot(c, c).real)) <= 1e-5
    ys = sample_indices(n, 23, 4096)
    got = qs.amplitudes(st, ys).astype(np.complex128)
    ref = closed.qft_wht_sparse(n, idx, c, closed.perm_source(n, perm, ys))
    assert rel_err(got, ref) <= REL["c64"], rel_err(got, ref)
    # index tags through the block alone
    t = st.tensor()
    chunk = 1 << 26
    for s in range(0, 1 << n, chunk):
        i = torch.arange(s, s + chunk, dtype=torch.int64, device="cuda")
        t[s:s + chunk] = torch.complex((i & ((1 << 24) - 1)).to(torch.float32), (i >> 24).to(torch.float32))
    qs.apply(st, qs.Plan(n, perm))
    ys = sample_indices(n, 29, 65536)
    src = closed.perm_source(n, perm, ys)
    want = ((src & np.uint64((1 << 24) - 1)).astype(np.float32)
            + 1j * (src >> np.uint64(24)).astype(np.float32)).astype(np.complex64)
    assert np.array_equal(qs.amplitudes(st, ys), want)
