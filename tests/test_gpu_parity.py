"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (floating point): state infidelity <= 1e-10 in complex64 and <= 1e-24
in complex128 (normalised, cancellation-free form), element-wise amplitude
agreement to a tolerance derived from float32 rounding; permutations are
bit-exact.  Inputs are seeded; the oracle starts from the device-rounded
input values.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed, metrics, statevec as sv

pytestmark = pytest.mark.gpu

INF64 = 1e-10
INF128 = 1e-24


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


def start(qs, n, dtype, seed=12):
    psi0 = W.gaussian_state(n, seed)
    nd = np.complex64 if dtype == "c64" else np.complex128
    psi0 = psi0.astype(nd)
    st = qs.State(n, dtype, init=None)
    st.upload(psi0)
    return st, psi0.astype(np.complex128)


def compare(qs, st, ref, dtype, n):
    got = st.download().astype(np.complex128)
    inf = metrics.infidelity(got, ref)
    bar = INF64 if dtype == "c64" else INF128
    assert inf <= bar, (n, dtype, inf)
    # element-wise: float32 rounding per operation, relative to the typical amplitude
    amp = 1.0 / math.sqrt(1 << n)
    atol = (5e-6 if dtype == "c64" else 1e-13) * amp * max(1.0, math.sqrt(n))
    assert np.max(np.abs(got - ref)) <= atol * 20, np.max(np.abs(got - ref)) / amp
    return inf


# ------------------------------------------------------------------ config 1: 12q QFT
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["plain", "fused"])
def test_qft12_gate_by_gate_and_fused(qs, dtype, mode):
    n = 12
    st, psi0 = start(qs, n, dtype)
    stream = W.qft_stream(n)
    if mode == "plain":
        qs.apply_gates(st, stream)
    else:
        qs.apply(st, qs.Plan(n, stream))
    ref = sv.run(psi0, n, stream)
    compare(qs, st, ref, dtype, n)
    assert abs(qs.norm2(st) - metrics.norm2(ref)) < (1e-6 if dtype == "c64" else 1e-14)


# ------------------------------------------------------------------ mixed streams
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (5, 4), (9, 5), (13, 6), (14, 7), (17, 8)])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_random_streams_plain_and_fused(qs, n, seed, dtype):
    kinds = None if n >= 2 else ("H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ", "P", "U")
    stream = W.random_stream(n, 150, seed, kinds)
    ref = None
    for mode in ("plain", "fused"):
        st, psi0 = start(qs, n, dtype, seed)
        if ref is None:
            ref = sv.run(psi0, n, stream)
        if mode == "plain":
            qs.apply_gates(st, stream)
        else:
            qs.apply(st, qs.Plan(n, stream))
        compare(qs, st, ref, dtype, n)


@pytest.mark.parametrize("tile_bits", [5, 8, 13, 14])
def test_tile_geometries(qs, tile_bits):
    n = 18
    stream = W.qft_stream(n) + W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 2, h_layer=False) + W.wht_stream(n)
    st, psi0 = start(qs, n, "c64", 3)
    plan = qs.Plan(n, stream, max_tile_bits=tile_bits)
    qs.apply(st, plan)
    compare(qs, st, sv.run(psi0, n, stream), "c64", n)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("case", ["approx2", "approx5", "adjacent", "adjacent_then_full"])
def test_approximate_and_register_qfts(qs, dtype, case):
    # stages whose bases differ (approximate QFT: stage p reads bits [p - d, p);
    # QFTs on neighbouring registers) share tile rounds; each computes its own
    # group twiddle
    n = 16
    if case.startswith("approx"):
        stream = W.qft_register_stream(range(n), int(case[-1]))
    else:
        hi, lo = W.qft_register_stream(range(7)), W.qft_register_stream(range(7, n))
        stream = lo + hi + (W.qft_stream(n) if case == "adjacent_then_full" else [])
    for tile_bits in (13, 7):
        st, psi0 = start(qs, n, dtype, 8)
        qs.apply(st, qs.Plan(n, stream, max_tile_bits=tile_bits))
        compare(qs, st, sv.run(psi0, n, stream), dtype, n)


def test_multi_qubit_and_controlled(qs):
    n = 11
    rng = np.random.default_rng(4)
    stream = (W.wht_stream(n) + [W.G("MCZ", 0, 3, 7), W.G("MCP", 1, 2, 9, 10, theta=0.3),
                                 W.G("UNITARY", 5, 1, 8, mat=W.random_unitary(8, rng)),
                                 W.G("UNITARY", 2, 6, mat=W.random_unitary(4, rng)),
                                 W.G("CU", 4, 0, mat=W.random_unitary(2, rng))] + W.random_stream(n, 40, 9))
    for mode in ("plain", "fused"):
        st, psi0 = start(qs, n, "c128", 5)
        if mode == "plain":
            qs.apply_gates(st, stream)
        else:
            qs.apply(st, qs.Plan(n, stream))
        compare(qs, st, sv.run(psi0, n, stream), "c128", n)


# ------------------------------------------------------------------ permutations (bit-exact)
@pytest.mark.parametrize("n", [2, 7, 12, 20])
def test_gf2_gather_bit_exact(qs, n):
    stream = W.random_perm_block(n, 200, 31)
    tag = W.index_tag_state(n).astype(np.complex64)
    for mode in ("plain", "fused"):
        st = qs.State(n, "c64", init=None)
        st.upload(tag)
        if mode == "plain":
            qs.apply_gates(st, stream)
        else:
            qs.apply(st, qs.Plan(n, stream))
        got = st.download()
        src = closed.perm_source(n, stream, np.arange(1 << n, dtype=np.uint64)).astype(np.int64)
        assert np.array_equal(got, tag[src]), mode


def test_ghz(qs):
    n = 16
    st = qs.State(n, "c64")
    qs.apply(st, qs.Plan(n, W.ghz_stream(n)))
    a = qs.amplitudes(st, [0, (1 << n) - 1, 1, 12345])
    assert np.allclose(a[:2], 1 / math.sqrt(2), atol=1e-7) and np.all(a[2:] == 0)


def test_grover_success(qs):
    n, k = 12, 8
    marked = 0b101100111010
    st = qs.State(n, "c128")
    qs.apply(st, qs.Plan(n, W.grover_stream(n, marked, k)))
    th = math.asin(1 / math.sqrt(1 << n))
    p = abs(qs.amplitudes(st, [marked])[0]) ** 2
    assert abs(p - math.sin((2 * k + 1) * th) ** 2) < 1e-12


# ------------------------------------------------------------------ reductions
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_expectations_norm_overlap(qs, dtype):
    n = 13
    st, psi = start(qs, n, dtype, 21)
    terms = W.xxz_terms(n, 0.5) + W.z_terms(n) + W.x_terms(n) + [(0.7, 0, 0), W.pauli(0.3, {0: "Y", 5: "X", 12: "Z"})]
    tot, per = qs.expect(st, terms, per_term=True)
    ref = sv.expect_terms(psi, n, terms)
    tol = 1e-7 if dtype == "c64" else 1e-13
    assert np.max(np.abs(per - ref)) < tol
    assert abs(tot - ref.sum()) < tol * len(terms)
    assert abs(qs.norm2(st) - metrics.norm2(psi)) < 1e-12
    st2, psi2 = start(qs, n, dtype, 22)
    ov = qs.overlap(st, st2)
    assert abs(ov - np.vdot(psi, psi2)) < 1e-12
    assert abs(qs.infidelity(st, st2) - metrics.infidelity(psi, psi2)) < 1e-12
    assert qs.infidelity(st, st) < 1e-28


def test_xxz_closed_forms_on_device(qs):
    n = 20
    terms = W.xxz_terms(n, 0.5)
    assert abs(qs.expect(qs.State(n, "c128"), terms) - 0.5 * (n - 1)) < 1e-12
    assert abs(qs.expect(qs.State(n, "c128", init="plus"), terms) - (n - 1)) < 1e-11
    neel = int("01" * (n // 2), 2)
    assert abs(qs.expect(qs.State(n, "c128").set_basis(neel), terms) + 0.5 * (n - 1)) < 1e-12


def test_reductions_are_deterministic(qs):
    n = 22
    st, _ = start(qs, n, "c64", 2)
    a = [qs.norm2(st) for _ in range(3)]
    b = [qs.expect(st, W.xxz_terms(n, 0.5)) for _ in range(3)]
    assert len(set(a)) == 1 and len(set(b)) == 1


# ------------------------------------------------------------------ invariants
def test_plan_then_inverse_returns_input(qs):
    n = 15
    stream = W.random_stream(n, 200, 13)
    st, psi0 = start(qs, n, "c128", 13)
    qs.apply(st, qs.Plan(n, stream))
    qs.apply(st, qs.Plan(n, sv.inverse_stream(stream)))
    assert metrics.infidelity(st.download(), psi0) < INF128


def test_error_paths_do_not_touch_the_state(qs):
    n = 6
    st, psi0 = start(qs, n, "c64", 1)
    with pytest.raises(qs.QsError):
        qs.apply(st, qs.Plan(7, W.wht_stream(7)))
    with pytest.raises(qs.QsError):
        qs.apply_gates(st, [W.G("H", 0), W.G("CNOT", 2, 2)])
    p = qs.Plan(n, [W.G("RX", 0, param=0)], n_params=1)
    with pytest.raises(qs.QsError):
        qs.apply(st, p)  # parameters not bound
    assert np.array_equal(st.download(), psi0.astype(np.complex64))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_empty_and_identity_plans(qs, dtype):
    """Degenerate plans: no gates, only identities, a gate and its inverse
    back to back; the state is returned unchanged (bit for bit where no
    arithmetic runs) and the fused norm falls back to a reduction."""
    n = 11
    st, psi0 = start(qs, n, dtype, 21)
    held = st.download().copy()
    for stream in ([], [W.G("I", q) for q in range(n)]):
        plan = qs.Plan(n, stream)
        assert plan.num_layers() == 0
        qs.apply(st, plan)
        qs.apply(st, plan.inverse())
        nrm = qs.apply_norm2(st, plan)
        assert np.array_equal(st.download(), held)
        h128 = held.astype(np.complex128)
        assert abs(nrm - float(np.vdot(h128, h128).real)) < 1e-12
    qs.apply(st, qs.Plan(n, [W.G("RX", 3, theta=0.4), W.G("RX", 3, theta=-0.4)]))
    tol = INF64 if dtype == "c64" else INF128
    assert metrics.infidelity(st.download(), held.astype(np.complex128)) <= tol


# ------------------------------------------------------------------ rotation layers
# Rotation rounds run in factored form when every |tan| <= 8 (one multiply-add
# per component, the cosines in the pass's store scale) and unfactored
# otherwise; both forms, negative cosines and the fused diagonal-then-rotation
# round are exercised, forward and through the inverse plan.
ROT_ANGLES = {
    "small": lambda q: 0.05 + 0.01 * q,
    "wide": lambda q: -2.5 + 0.4 * q,
    "near_pi": lambda q: math.pi - 0.01 * (q + 1),
    "mixed": lambda q: [0.3, math.pi - 0.02, -1.1, 2.9, 0.7][q % 5],
}


@pytest.mark.parametrize("kind", ["RX", "RY"])
@pytest.mark.parametrize("angles", sorted(ROT_ANGLES))
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_rotation_layers_factored_and_plain_forms(qs, kind, angles, dtype):
    n = 16
    f = ROT_ANGLES[angles]
    stream = []
    for layer in range(3):
        stream += [W.G(kind, q, theta=f(q) * (1.0 + 0.1 * layer)) for q in range(n)]
        stream += [W.G("RZZ", q, q + 1, theta=0.3 + 0.05 * layer) for q in range(n - 1)]
    stream += [W.G(kind, q, theta=f(n - 1 - q)) for q in range(n)]
    st, psi0 = start(qs, n, dtype)
    plan = qs.Plan(n, stream, max_tile_bits=8)
    qs.apply(st, plan)
    ref = sv.run(psi0, n, stream)
    compare(qs, st, ref, dtype, n)
    assert abs(qs.norm2(st) - metrics.norm2(ref)) < (1e-6 if dtype == "c64" else 1e-13)
    qs.apply(st, plan.inverse())
    compare(qs, st, psi0, dtype, n)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("dl,bal", [(0, 0), (-1, 0), (-1, -1), (4, 0)])
def test_tfim_diagonal_pass_options_match_oracle(qs, dtype, dl, bal):
    n = 18
    stream = W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 6)
    st, psi0 = start(qs, n, dtype)
    qs.apply(st, qs.Plan(n, stream, max_tile_bits=10, diag_low_bits=dl, balance_passes=bal))
    compare(qs, st, sv.run(psi0, n, stream), dtype, n)


def test_long_rotation_runs_keep_the_norm(qs):
    # 60 Strang steps at 20 qubits in complex64: the factored rotations' scales
    # are rounded with the running norm compensation
    n = 20
    stream = W.tfim_strang_stream(n, 1.0, 0.9, 0.07, 60)
    st, _ = start(qs, n, "c64")
    before = qs.norm2(st)
    qs.apply(st, qs.Plan(n, stream))
    assert abs(qs.norm2(st) / before - 1.0) < 2e-6


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_single_qubit_round_factorisations(qs, dtype):
    """Layers of single-qubit gates whose fused 2x2 matrices sit at the edges
    of the tile rounds' D2 [[1, -t], [t, 1]] D1 form: pure phases (t = 0),
    X-like matrices (no factorisation: the plain matrix round), |t| just below
    and above the factored bound 8, Hadamards (scaled unitaries), RY near pi,
    RY then RZ (D1 all ones), RZ then RY (D2 all ones) and Haar unitaries
    (both tables), three layers deep, against the oracle."""
    n = 14
    rng = np.random.default_rng(21)
    t8 = 2.0 * math.atan(8.0)
    per_qubit = [
        [W.G("RZ", 0, theta=0.7), W.G("S", 0), W.G("T", 0)],
        [W.G("X", 0), W.G("RZ", 0, theta=0.3)],
        [W.G("RY", 0, theta=t8 - 1e-3)],
        [W.G("RY", 0, theta=t8 + 1e-3)],
        [W.G("H", 0)],
        [W.G("RY", 0, theta=math.pi - 1e-4), W.G("RZ", 0, theta=-1.1)],
        [W.G("RY", 0, theta=0.4), W.G("RZ", 0, theta=1.3)],
        [W.G("RZ", 0, theta=-0.6), W.G("RY", 0, theta=2.2)],
        [W.G("U", 0, mat=W.random_unitary(2, rng))],
        [W.G("SX", 0), W.G("P", 0, theta=0.9)],
        [W.G("Y", 0)],
        [W.G("RX", 0, theta=1.7), W.G("RZ", 0, theta=0.2)],
        [W.G("U", 0, mat=W.random_unitary(2, rng)), W.G("H", 0)],
        [W.G("RY", 0, theta=-2.9)],
    ]
    stream = []
    for layer in range(3):
        for q in range(n):
            for g in per_qubit[(q + 5 * layer) % len(per_qubit)]:
                mat = None if g.mat is None else np.array(g.mat).reshape(2, 2)
                stream.append(W.G(g.name, q, theta=g.theta, mat=mat))
        stream.append(W.G("CNOT", layer, layer + 7))
    st, psi0 = start(qs, n, dtype, 4)
    plan = qs.Plan(n, stream, window_k=-1)  # structured tile rounds, no dense windows
    assert all(l["kind"] != "dense" for l in plan.describe()["layers"])
    qs.apply(st, plan)
    compare(qs, st, sv.run(psi0, n, stream), dtype, n)
